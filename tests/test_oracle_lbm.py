"""Pins of the oracle's lattice Boltzmann part (Section 2.1, eqs 5-11).

Each check is fixed by the mathematics, not by re-running the oracle's own
formula: moments of the equilibrium (eq 6), the mass and momentum budget of
the Guo forcing scheme (eqs 5, 7, 11), uniform flow, the analytic
body-force Poiseuille profile with halfway bounce-back walls, and the
viscous decay rate of a shear wave (the viscosity-relaxation relation).
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

# eq 8
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def sim(nx, ny, bc=W.FULLY_PERIODIC, tau=0.8, G=(0.0, 0.0), inflow=(0.0, 0.0), init=(1.0, 0.0, 0.0)):
    return OracleSim(nx, ny, bc, tau, W.COS4, 2.6, G, inflow, init)


def moment(f, a, b):
    return np.einsum("q,q,qij->ij", a, b, f)


def test_equilibrium_moments(oracle_lib):
    rng = np.random.default_rng(0)
    nx, ny = 11, 7
    rho = 1 + 0.05 * rng.standard_normal((ny, nx))
    ux = 0.05 * rng.standard_normal((ny, nx))
    uy = 0.05 * rng.standard_normal((ny, nx))
    s = sim(nx, ny)
    s.init_equilibrium(ux, uy, rho)
    f = s.populations()
    one = np.ones(9)
    assert np.allclose(moment(f, one, one), rho, rtol=0, atol=1e-15)
    assert np.allclose(moment(f, EX, one), rho * ux, rtol=0, atol=1e-16)
    assert np.allclose(moment(f, EY, one), rho * uy, rtol=0, atol=1e-16)
    # second moments: rho (u u + I/3)
    assert np.allclose(moment(f, EX, EX), rho * (ux * ux + 1 / 3), rtol=0, atol=1e-15)
    assert np.allclose(moment(f, EX, EY), rho * ux * uy, rtol=0, atol=1e-16)
    assert np.allclose(moment(f, EY, EY), rho * (uy * uy + 1 / 3), rtol=0, atol=1e-15)


def test_mass_and_momentum_budget_with_body_force(oracle_lib):
    # Guo scheme: per node, sum_q A' = rho and sum_q e_q A' = m + f (so the
    # total momentum grows by exactly N G per step on a periodic grid)
    rng = np.random.default_rng(1)
    nx, ny = 23, 17
    G = (3e-5, -2e-5)
    s = sim(nx, ny, G=G, tau=0.63)
    ux = 0.04 * np.sin(2 * np.pi * np.arange(ny) / ny)[:, None] * np.ones((1, nx))
    uy = 0.02 * rng.standard_normal((ny, nx))
    rho = 1 + 0.01 * rng.standard_normal((ny, nx))
    s.init_equilibrium(ux, uy, rho)
    one = np.ones(9)
    for _ in range(5):
        r, us, vs = s.macroscopic()         # moments of the streamed populations
        mx = r * us - 0.5 * G[0]
        my = r * vs - 0.5 * G[1]
        f0 = s.populations()
        s.step(1)
        f1 = s.populations()
        assert np.allclose(moment(f1, one, one), r, rtol=0, atol=2e-15)
        assert np.allclose(moment(f1, EX, one), mx + G[0], rtol=0, atol=2e-16)
        assert np.allclose(moment(f1, EY, one), my + G[1], rtol=0, atol=2e-16)
        assert abs(f1.sum() - f0.sum()) < 1e-12
        px0, px1 = moment(f0, EX, one).sum(), moment(f1, EX, one).sum()
        assert abs(px1 - px0 - nx * ny * G[0]) < 1e-13


@pytest.mark.parametrize("bc", [W.FULLY_PERIODIC, W.CHANNEL])
def test_uniform_flow_stays_uniform(oracle_lib, bc):
    u0 = (0.03, 0.0) if bc == W.CHANNEL else (0.03, -0.01)
    s = sim(40, 20, bc=bc, inflow=u0, init=(1.0,) + u0)
    f0 = s.populations()
    s.step(50)
    assert np.max(np.abs(s.populations() - f0)) < 1e-15


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.5, 0.5 + np.sqrt(3) / 4])
def test_poiseuille_bounce_back(oracle_lib, tau):
    # walls at y = -1/2 and y = H - 1/2 (halfway bounce-back); with y = j + 1/2
    # the steady discrete solution is u = G/(2 nu) y (H - y) + G (16 tau^2 - 16 tau + 1)/(24 nu)
    H, G = 16, 1e-6
    nu = (tau - 0.5) / 3
    s = sim(4, H, bc=(W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), tau=tau, G=(G, 0.0))
    steps = int(40 * H * H / (np.pi ** 2 * nu)) + 1000
    s.step(steps)
    _, u, v = s.macroscopic()
    y = np.arange(H) + 0.5
    exact = G / (2 * nu) * y * (H - y) + G * (16 * tau * tau - 16 * tau + 1) / (24 * nu)
    # u* includes G/2; the collision velocity is u* (no IB force here), so compare u*
    assert np.max(np.abs(u[:, 1] - exact)) < 1e-9 * np.max(exact)
    assert np.max(np.abs(v)) < 1e-10 * np.max(exact)
    # curvature -G/nu exactly
    d2 = u[2:, 1] - 2 * u[1:-1, 1] + u[:-2, 1]
    assert np.allclose(d2, -G / nu, rtol=1e-8, atol=0)


def test_shear_wave_viscosity(oracle_lib):
    # u_x = A sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3
    ny, tau = 64, 0.8
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / ny
    s = sim(4, ny, tau=tau)
    y = np.arange(ny)
    ux = 1e-3 * np.sin(k * y)[:, None] * np.ones((1, 4))
    s.init_equilibrium(ux, np.zeros_like(ux))

    def amp():
        _, u, _ = s.macroscopic()
        return 2 * np.mean(u[:, 0] * np.sin(k * y))

    s.step(200)
    a0 = amp()
    s.step(2000)
    a1 = amp()
    rate = -np.log(a1 / a0) / 2000
    assert abs(rate / (nu * k * k) - 1) < 2e-3
