"""The oracle's rigid body motion (eq 4 for a rigid body: the surface
moves with the fluid it carries, U_l = V + omega x (X_l - c)).

Pins: the closed-form kinematics after n steps; a body carried along by a
uniform flow at the flow's own velocity feels no force and leaves the flow
exactly as it was; a body set in motion with zero velocity is a fixed body;
the fluid's momentum changes each step by exactly minus the force on the
bodies (eq 27), with bodies translating and turning.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])[:, None, None]
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])[:, None, None]


def test_closed_form_kinematics():
    o = OracleSim(64, 64, W.FULLY_PERIODIC, 0.8, W.ROMA3, 1.9)
    b = W.cylinder_body(30.2, 29.7, 10.0, 31)
    o.add_body(b.xy, None, b.cx, b.cy, b.ds)
    V, om = (0.013, -0.007), 0.004
    o.set_body_motion(0, V[0], V[1], om)
    n = 37
    o.step(n)
    st = o.body_state(0)
    c = np.array([b.cx + n * V[0], b.cy + n * V[1]])
    assert np.max(np.abs(st[:2] - c)) < 1e-12 and abs(st[2] - n * om) < 1e-14
    r = b.xy - [b.cx, b.cy]
    R = np.array([[np.cos(n * om), -np.sin(n * om)], [np.sin(n * om), np.cos(n * om)]])
    assert np.max(np.abs(o.marker_positions() - (c + r @ R.T))) < 1e-12


def test_marker_velocity_is_the_rigid_field():
    """Read back through the force of a comoving uniform flow: U_l must be
    V + omega x (X_l - c); checked on the interpolated direct force."""
    o = OracleSim(64, 64, W.FULLY_PERIODIC, 0.8, W.ROMA3, 1.9, init=(1.0, 0.0, 0.0))
    b = W.cylinder_body(30.2, 29.7, 10.0, 31)
    o.add_body(b.xy, None, b.cx, b.cy, b.ds)
    om = 0.003
    o.set_body_motion(0, 0.0, 0.0, om)
    o.step(1)
    md = o.marker_data()  # fluid at rest: F_l = 2 rho_l U_l
    xy0 = b.xy - [b.cx, b.cy]
    U = np.stack([-om * xy0[:, 1], om * xy0[:, 0]], axis=1)
    assert np.max(np.abs(md["Fx"] - 2 * md["rho"] * U[:, 0])) < 1e-15
    assert np.max(np.abs(md["Fy"] - 2 * md["rho"] * U[:, 1])) < 1e-15


@pytest.mark.parametrize("kind", [W.ROMA3, W.COS4])
def test_a_body_carried_by_a_uniform_flow_feels_nothing(kind):
    V = (0.031, -0.012)
    o = OracleSim(64, 48, W.FULLY_PERIODIC, 0.8, kind, 1.9, init=(1.0, *V))
    b = W.cylinder_body(20.3, 22.6, 9.0, 28)
    o.add_body(b.xy, None, b.cx, b.cy, b.ds)
    o.set_body_motion(0, *V, 0.0)
    f0 = o.populations()
    for _ in range(60):
        o.step(1)
        assert np.max(np.abs(o.forces())) < 1e-13
    assert np.max(np.abs(o.populations() - f0)) < 1e-13
    assert abs(o.body_state(0)[0] - (20.3 + 60 * V[0])) < 1e-12


def test_zero_motion_is_a_fixed_body():
    c = W.random_case(60, nx=60, ny=50, kind=W.PESKIN4, bc=W.FULLY_PERIODIC, n_bodies=2, moving=False)
    runs = []
    for move in (False, True):
        o = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
        for b in c.bodies:
            o.add_body(b.xy, None, b.cx, b.cy, b.ds)
        if move:
            o.set_body_motion(1, 0.0, 0.0, 0.0)
        o.step(10)
        runs.append(o.populations())
    assert np.max(np.abs(runs[0] - runs[1])) < 1e-14


@pytest.mark.parametrize("bc", [W.FULLY_PERIODIC, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL)])
def test_fluid_momentum_balances_the_body_forces(bc):
    """Guo forcing adds the spread force to the fluid's momentum and the
    force on the bodies is minus that force (eq 27): with no body force and
    a fully periodic grid the x-momentum changes by -sum F_x each step.
    Mass is conserved with walls too."""
    o = OracleSim(72, 56, bc, 0.75, W.ROMA3, 1.9, init=(1.0, 0.0, 0.0))
    b1 = W.cylinder_body(25.3, 27.1, 10.0, 31)
    b2 = W.cylinder_body(50.1, 30.4, 8.0, 25)
    o.add_body(b1.xy, None, b1.cx, b1.cy, b1.ds)
    o.add_body(b2.xy, None, b2.cx, b2.cy, b2.ds)
    o.set_body_motion(0, 0.02, 0.004, 0.002)
    o.set_body_motion(1, -0.01, 0.0, -0.003)
    f = o.populations()
    for _ in range(20):
        px, mass = (EX * f).sum(), f.sum()
        o.step(1)
        f = o.populations()
        F = o.forces()
        assert abs(f.sum() - mass) < 1e-12
        if bc == W.FULLY_PERIODIC:
            assert abs((EX * f).sum() - px + F[:, 0].sum()) < 1e-12
