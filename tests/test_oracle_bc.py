"""The oracle's far-field boundaries of the cylinder runs (Section 5.2).

Free-slip walls (du_x/dy = 0, u_y = 0 at the top and bottom) are realised as
a specular reflection halfway between the edge row and the wall; the
convective outlet advects the ghost column with the inflow speed U,
implicit upwind: phi_N(t+1) = (phi_N(t) + U phi_{N-1}(t+1)) / (1 + U).
Neither realisation is printed in the paper; the pins below fix them by
what the continuous conditions imply:

* method of images: a free-slip channel of height ny evolves exactly as the
  lower half of a periodic channel of height 2 ny holding the mirror-image
  flow (and the mirror-image bodies);
* closed forms: uniform flow along free-slip walls is a fixed point, and a
  uniform body force accelerates the whole channel uniformly, u = (n + 1/2) G;
* conservation: mass and x-momentum, exactly, with no body force;
* the convective outlet: a uniform inflow is a fixed point; with U = 0 the
  ghost column is frozen; d(ghost)/dU at U = 0 equals the difference of the
  new column nx-2 and the old ghost (the discrete equation's first-order
  term); steady states equal those of the zero-gradient outlet.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

SLIP_Y = (W.PERIODIC, W.PERIODIC, W.FREE_SLIP_WALL, W.FREE_SLIP_WALL)
MIRROR = [0, 1, 4, 3, 2, 8, 7, 6, 5]  # q -> the direction with (e_x, -e_y), D2Q9 order of eq 8


def random_fields(rng, nx, ny, amp=0.02):
    rho = 1.0 + 0.5 * amp * rng.uniform(-1, 1, size=(ny, nx))
    ux = amp * rng.uniform(-1, 1, size=(ny, nx))
    uy = amp * rng.uniform(-1, 1, size=(ny, nx))
    return rho, ux, uy


@pytest.mark.parametrize("kind", [W.ROMA3, W.COS4])
def test_free_slip_is_the_mirror_image_of_a_periodic_channel(kind):
    nx, ny, n = 24, 14, 30
    rng = np.random.default_rng(3)
    rho, ux, uy = random_fields(rng, nx, ny)
    G = (2e-5, 0.0)
    body = W.cylinder_body(10.3, 6.2, 5.0, n=13)
    uv = rng.uniform(-0.01, 0.01, size=(13, 2))

    s = OracleSim(nx, ny, SLIP_Y, 0.8, kind, 1.9, G)
    s.add_body(body.xy, uv, body.cx, body.cy, body.ds)
    s.init_equilibrium(ux, uy, rho)

    d = OracleSim(nx, 2 * ny, W.FULLY_PERIODIC, 0.8, kind, 1.9, G)
    d.add_body(body.xy, uv, body.cx, body.cy, body.ds)
    mxy = np.stack([body.xy[:, 0], (2 * ny - 1) - body.xy[:, 1]], axis=1)
    muv = np.stack([uv[:, 0], -uv[:, 1]], axis=1)
    d.add_body(mxy, muv, body.cx, (2 * ny - 1) - body.cy, body.ds)
    d.init_equilibrium(np.vstack([ux, ux[::-1]]), np.vstack([uy, -uy[::-1]]), np.vstack([rho, rho[::-1]]))

    for step in range(n):
        s.step(1)
        d.step(1)
        fs, fd = s.populations(), d.populations()
        assert np.max(np.abs(fd[:, :ny] - fs)) < 1e-14, step
        # the upper half stays the mirror image
        assert np.max(np.abs(fd[MIRROR, ny:][:, ::-1] - fs)) < 1e-14, step
    Fs, Fd = s.forces(), d.forces()
    assert np.max(np.abs(Fd[0] - Fs[0])) < 1e-12 * np.max(np.abs(Fs))
    assert np.max(np.abs(Fd[1] * [1, -1, -1] - Fs[0])) < 1e-12 * np.max(np.abs(Fs))


def test_uniform_flow_along_free_slip_walls_is_a_fixed_point():
    nx, ny = 20, 10
    for bc, fixed in ((SLIP_Y, True), ((W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), False)):
        s = OracleSim(nx, ny, bc, 0.7, W.ROMA3, 1.9, init=(1.0, 0.05, 0.0))
        f0 = s.populations()
        s.step(200)
        moved = np.max(np.abs(s.populations() - f0))
        assert (moved < 1e-15) == fixed, (bc, moved)


def test_body_force_accelerates_a_free_slip_channel_uniformly():
    """Guo forcing adds G to the momentum of every node each step; with
    free-slip walls nothing opposes it, so u = (n + 1/2) G / rho everywhere."""
    nx, ny, G = 16, 12, 3e-6
    s = OracleSim(nx, ny, SLIP_Y, 0.9, W.ROMA3, 1.9, (G, 0.0))
    for n in (1, 10, 100):
        s.step(n - s.steps)
        rho, ux, uy = s.macroscopic()
        assert np.max(np.abs(rho - 1.0)) < 1e-13
        assert np.max(np.abs(ux - (n + 0.5) * G)) < 1e-13
        assert np.max(np.abs(uy)) < 1e-14


def test_free_slip_conserves_mass_and_x_momentum():
    nx, ny = 30, 16
    rng = np.random.default_rng(4)
    rho, ux, uy = random_fields(rng, nx, ny, amp=0.03)
    s = OracleSim(nx, ny, SLIP_Y, 0.75, W.ROMA3, 1.9)
    s.init_equilibrium(ux, uy, rho)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])[:, None, None]
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])[:, None, None]
    f = s.populations()
    m0, px0, py0 = f.sum(), (ex * f).sum(), (ey * f).sum()
    drift_y = 0.0
    for _ in range(40):
        s.step(1)
        f = s.populations()
        assert abs(f.sum() - m0) < 1e-14 * m0
        assert abs((ex * f).sum() - px0) < 1e-14 * m0
        drift_y = max(drift_y, abs((ey * f).sum() - py0))
    assert drift_y > 1e-6  # the walls do exchange y-momentum


def far_field(nx, ny, U, tau=0.8, G=(0.0, 0.0), outlet=W.CONVECTIVE_OUTLET):
    return OracleSim(nx, ny, (W.VELOCITY_INLET, outlet, W.FREE_SLIP_WALL, W.FREE_SLIP_WALL), tau, W.ROMA3,
                     1.9, G, (U, 0.0), (1.0, U, 0.0))


def test_uniform_inflow_is_a_fixed_point_of_the_far_field_boundaries():
    s = far_field(30, 12, 0.05)
    f0 = s.populations()
    s.step(300)
    assert np.max(np.abs(s.populations() - f0)) < 1e-15


def test_convective_outlet_ghost_is_frozen_at_zero_speed():
    nx, ny = 24, 10
    rng = np.random.default_rng(5)
    rho, ux, uy = random_fields(rng, nx, ny)
    s = far_field(nx, ny, 0.0)
    s.init_equilibrium(ux, uy, rho)
    g0 = s.populations()[:, :, -1].copy()
    s.step(25)
    f = s.populations()
    assert np.array_equal(f[:, :, -1], g0)
    assert np.max(np.abs(f[:, :, -2] - g0)) > 1e-4


def test_convective_outlet_first_order_in_the_speed():
    """phi_N(t+1) - phi_N(t) = U (phi_{N-1}(t+1) - phi_N(t)) + O(U^2)."""
    nx, ny = 24, 10
    rng = np.random.default_rng(6)
    rho, ux, uy = random_fields(rng, nx, ny)
    out = {}
    for U in (0.0, 1e-6, 2e-6):
        s = far_field(nx, ny, U)
        s.init_equilibrium(ux, uy, rho)
        old = s.populations()[:, :, -1].copy()
        s.step(1)
        f = s.populations()
        out[U] = (f[:, :, -1], f[:, :, -2])
    # column nx-2 does not see the inflow speed after one step
    assert np.array_equal(out[0.0][1], out[1e-6][1])
    expect = out[0.0][1] - old
    for U in (1e-6, 2e-6):
        deriv = (out[U][0] - out[0.0][0]) / U   # = expect / (1 + U) exactly
        assert np.max(np.abs(deriv - expect)) < 2 * U * np.max(np.abs(expect)) + 1e-9


def test_convective_and_zero_gradient_outlets_share_steady_states():
    nx, ny, U = 48, 20, 0.04
    body = W.cylinder_body(14.3, 10.2, 6.0)
    runs = []
    for outlet in (W.CONVECTIVE_OUTLET, W.ZERO_GRADIENT_OUTLET):
        s = far_field(nx, ny, U, tau=0.9, outlet=outlet)
        s.add_body(body.xy, None, body.cx, body.cy, body.ds)
        s.step(6000)
        a = s.populations()
        s.step(1)
        b = s.populations()
        assert np.max(np.abs(b - a)) < 1e-13, outlet   # steady
        runs.append(b)
    # at a steady state the convective ghost equals column nx-2
    assert np.max(np.abs(runs[0][:, :, -1] - runs[0][:, :, -2])) < 1e-12
    # so the steady equations are those of the zero-gradient outlet; they
    # leave the mean density free (f -> c f maps steady states to steady
    # states: the collision, the direct force 2 rho (U - u) and both ghost
    # columns are homogeneous of degree one), so the two runs agree up to c
    c = runs[0][:, :, 1:-1].sum() / runs[1][:, :, 1:-1].sum()
    assert abs(c - 1.0) > 1e-4
    assert np.max(np.abs(runs[0] - c * runs[1])) < 1e-12
